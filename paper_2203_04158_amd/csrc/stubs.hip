// Entry points whose implementation has not landed yet report EUNSUPPORTED.
#include "common.hpp"

struct LearnedModel {};

void learned_free(LearnedModel *m) { delete m; }
uint64_t learned_bytes(const LearnedModel *) { return 0; }

mbr_status rank_learned_launch(const mbr_ranker *, const void *, uint64_t, uint32_t *, hipStream_t) {
    MBR_FAIL(MBR_EUNSUPPORTED, "learned ranking not built");
}

extern "C" {
mbr_status mbr_learned_train(const mbr_sector *, const mbr_learned_opts *, const mbr_ranker *,
                             mbr_ranker **, void *) {
    MBR_FAIL(MBR_EUNSUPPORTED, "learned index not built");
}
mbr_status mbr_learned_max_error(const mbr_ranker *, uint64_t *, int32_t *) {
    MBR_FAIL(MBR_EUNSUPPORTED, "learned index not built");
}
mbr_status mbr_learned_params(const mbr_ranker *, float *, void *) {
    MBR_FAIL(MBR_EUNSUPPORTED, "learned index not built");
}
mbr_status mbr_mlp_forward(const float *, const uint32_t *, int32_t, float *, void *) {
    MBR_FAIL(MBR_EUNSUPPORTED, "learned index not built");
}
mbr_status mbr_mlp_gradients(const float *, const uint32_t *, const float *, int32_t, float *,
                             float *, void *) {
    MBR_FAIL(MBR_EUNSUPPORTED, "learned index not built");
}
}
