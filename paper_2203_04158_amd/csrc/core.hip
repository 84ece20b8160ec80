// Error reporting, binomial tables, handle bookkeeping and the rank dispatcher.
#include <cstdarg>
#include <mutex>

#include "common.hpp"

namespace mbr {

static thread_local std::string g_err;

void set_error(const char *fmt, ...) {
    char buf[1024];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    g_err = buf;
}

void clear_error() { g_err.clear(); }

mbr_status upload(DevBuf &b, const void *host, size_t bytes, hipStream_t stream) {
    MBR_TRY(b.alloc(bytes));
    if (bytes) {
        MBR_HIP(hipMemcpyAsync(b.p, host, bytes, hipMemcpyHostToDevice, stream));
        MBR_HIP(hipStreamSynchronize(stream));
    }
    return MBR_OK;
}

static uint64_t g_binom[65][65];
static std::once_flag g_binom_once;

static void binom_fill() {
    for (int n = 0; n <= 64; ++n) {
        g_binom[n][0] = 1;
        for (int k = 1; k <= 64; ++k)
            g_binom[n][k] = n == 0 ? 0 : g_binom[n - 1][k - 1] + g_binom[n - 1][k];
    }
}

uint64_t binom(int n, int k) {
    std::call_once(g_binom_once, binom_fill);
    if (n < 0 || k < 0 || n > 64 || k > 64) return 0;
    return g_binom[n][k];
}

static std::mutex g_dev_mutex;
static void *g_dev_binom[64] = {nullptr};

mbr_status device_binom(const uint64_t **d_table) {
    int dev = 0;
    MBR_HIP(hipGetDevice(&dev));
    if (dev < 0 || dev >= 64) MBR_FAIL(MBR_EUNSUPPORTED, "device index %d", dev);
    std::lock_guard<std::mutex> lk(g_dev_mutex);
    if (!g_dev_binom[dev]) {
        binom(0, 0);
        void *p = nullptr;
        MBR_HIP(hipMalloc(&p, sizeof g_binom));
        MBR_HIP(hipMemcpy(p, g_binom, sizeof g_binom, hipMemcpyHostToDevice));
        g_dev_binom[dev] = p;
    }
    *d_table = static_cast<const uint64_t *>(g_dev_binom[dev]);
    return MBR_OK;
}

int device_cu_count() {
    int dev = 0, cus = 0;
    if (hipGetDevice(&dev) != hipSuccess) return 256;
    if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess ||
        cus <= 0)
        return 256;
    return cus;
}

}  // namespace mbr

mbr_ranker::~mbr_ranker() {
    if (trie) trie_free(trie);
    if (btrie) bitmap_trie_free(btrie);
    if (learned) learned_free(learned);
}

extern "C" {

const char *mbr_status_str(mbr_status s) {
    switch (s) {
        case MBR_OK: return "ok";
        case MBR_EINVAL: return "invalid argument";
        case MBR_ENOMEM: return "out of memory";
        case MBR_EHIP: return "HIP runtime error";
        case MBR_ENOTSORTED: return "state list not sorted";
        case MBR_EDUP: return "state list has duplicates";
        case MBR_ERANGE: return "index or size out of range";
        case MBR_EUNSUPPORTED: return "unsupported";
        default: return "unknown status";
    }
}

const char *mbr_last_error(void) { return mbr::g_err.c_str(); }

int32_t mbr_version(void) { return 10100; }

mbr_status mbr_trie_bytes(const mbr_ranker *r, uint64_t *bytes) {
    if (!r || !bytes) MBR_FAIL(MBR_EINVAL, "null ranker or output");
    if (r->kind == MBR_RANKER_TRIE) *bytes = trie_bytes(r->trie);
    else if (r->kind == MBR_RANKER_BITMAP_TRIE) *bytes = r->btrie ? r->btrie->table.bytes : 0;
    else MBR_FAIL(MBR_EINVAL, "not a trie ranker (kind %d)", r->kind);
    return MBR_OK;
}

mbr_status mbr_ranker_info_get(const mbr_ranker *r, mbr_ranker_info *info) {
    if (!r || !info) MBR_FAIL(MBR_EINVAL, "null ranker or info");
    mbr_ranker_info o{};
    o.kind = r->kind;
    o.M = r->M;
    o.k = r->k;
    o.width_bits = r->width_bits;
    o.n_states = r->n_states;
    switch (r->kind) {
        case MBR_RANKER_STAGGERED:
        case MBR_RANKER_SPIN:
            o.bytes = r->stag.table.bytes;
            o.levels = r->stag.nch;
            break;
        case MBR_RANKER_TRIE:
            o.bytes = trie_bytes(r->trie);
            o.levels = trie_levels(r->trie);
            break;
        case MBR_RANKER_LEARNED:
            o.bytes = learned_bytes(r->learned);
            o.levels = 0;
            break;
        case MBR_RANKER_BITMAP_TRIE:
            o.bytes = r->btrie ? r->btrie->table.bytes : 0;
            o.levels = r->btrie ? r->btrie->H : 0;
            break;
        case MBR_RANKER_SAMPLED:
            o.bytes = learned_bytes(r->learned);
            o.levels = learned_levels(r->learned);
            break;
        case MBR_RANKER_BISECT:
            o.bytes = r->sector ? r->sector->states.bytes : 0;
            o.levels = 0;
            break;
        case MBR_RANKER_CNS:
            o.bytes = r->stag.table.bytes;
            o.levels = r->N;
            break;
        default: break;
    }
    *info = o;
    return MBR_OK;
}

mbr_status mbr_rank_batch(const mbr_ranker *r, const void *d_q, uint64_t n, uint32_t *d_rank,
                          void *stream) {
    if (!r) MBR_FAIL(MBR_EINVAL, "null ranker");
    if (n == 0) return MBR_OK;
    if (!d_q || !d_rank) MBR_FAIL(MBR_EINVAL, "null query or output pointer");
    if (n > (uint64_t)1 << 40) MBR_FAIL(MBR_ERANGE, "batch of %llu queries", (unsigned long long)n);
    hipStream_t s = mbr::as_stream(stream);
    switch (r->kind) {
        case MBR_RANKER_STAGGERED: return rank_staggered_launch(r, d_q, n, d_rank, s);
        case MBR_RANKER_SPIN: return rank_spin_launch(r, d_q, n, d_rank, s);
        case MBR_RANKER_TRIE: return rank_trie_launch(r, d_q, n, d_rank, s);
        case MBR_RANKER_BITMAP_TRIE: return rank_bitmap_trie_launch(r, d_q, n, d_rank, s);
        case MBR_RANKER_LEARNED:
        case MBR_RANKER_SAMPLED: return rank_learned_launch(r, d_q, n, d_rank, s);
        case MBR_RANKER_BISECT: return rank_bisect_launch(r, d_q, n, d_rank, s);
        case MBR_RANKER_CNS: return rank_cns_launch(r, d_q, n, d_rank, s);
        default: MBR_FAIL(MBR_EINVAL, "unknown ranker kind %d", r->kind);
    }
}

mbr_status mbr_rank_batch64(const mbr_ranker *r, const void *d_q, uint64_t n, uint64_t *d_rank,
                            void *stream) {
    if (!r) MBR_FAIL(MBR_EINVAL, "null ranker");
    if (n == 0) return MBR_OK;
    if (!d_q || !d_rank) MBR_FAIL(MBR_EINVAL, "null query or output pointer");
    if (n > (uint64_t)1 << 40) MBR_FAIL(MBR_ERANGE, "batch of %llu queries", (unsigned long long)n);
    if (r->kind != MBR_RANKER_STAGGERED)
        MBR_FAIL(MBR_EUNSUPPORTED, "64-bit ranks come from staggered rankers only");
    return rank_staggered_launch64(r, d_q, n, d_rank, mbr::as_stream(stream));
}

mbr_status mbr_ranker_destroy(mbr_ranker *r) {
    delete r;
    return MBR_OK;
}

}  // extern "C"
