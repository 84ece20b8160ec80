// Entry points whose implementation has not landed yet report EUNSUPPORTED.
#include "common.hpp"

struct TrieLevels {};
struct LearnedModel {};

void trie_free(TrieLevels *t) { delete t; }
uint64_t trie_bytes(const TrieLevels *) { return 0; }
int32_t trie_levels(const TrieLevels *) { return 0; }
void learned_free(LearnedModel *m) { delete m; }
uint64_t learned_bytes(const LearnedModel *) { return 0; }

mbr_status rank_trie_launch(const mbr_ranker *, const void *, uint64_t, uint32_t *, hipStream_t) {
    MBR_FAIL(MBR_EUNSUPPORTED, "trie ranking not built");
}
mbr_status rank_learned_launch(const mbr_ranker *, const void *, uint64_t, uint32_t *, hipStream_t) {
    MBR_FAIL(MBR_EUNSUPPORTED, "learned ranking not built");
}

extern "C" {
mbr_status mbr_build_trie(const mbr_sector *, int32_t, mbr_ranker **, void *) {
    MBR_FAIL(MBR_EUNSUPPORTED, "trie not built");
}
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
mbr_status mbr_hubbard_create(const mbr_hubbard_desc *, mbr_hubbard **, void *) {
    MBR_FAIL(MBR_EUNSUPPORTED, "not built");
}
mbr_status mbr_hubbard_dim(const mbr_hubbard *, uint64_t *, uint64_t *) { MBR_FAIL(MBR_EUNSUPPORTED, "not built"); }
mbr_status mbr_hubbard_apply(const mbr_hubbard *, const void *, void *, void *) { MBR_FAIL(MBR_EUNSUPPORTED, "not built"); }
mbr_status mbr_hubbard_destroy(mbr_hubbard *) { return MBR_OK; }
mbr_status mbr_lanczos_create(const mbr_hubbard *, const mbr_lanczos_opts *, mbr_lanczos **) { MBR_FAIL(MBR_EUNSUPPORTED, "not built"); }
mbr_status mbr_lanczos_start(mbr_lanczos *, const double *, void *) { MBR_FAIL(MBR_EUNSUPPORTED, "not built"); }
mbr_status mbr_lanczos_step(mbr_lanczos *, int32_t, void *) { MBR_FAIL(MBR_EUNSUPPORTED, "not built"); }
mbr_status mbr_lanczos_result(mbr_lanczos *, double *, int32_t *, void *) { MBR_FAIL(MBR_EUNSUPPORTED, "not built"); }
mbr_status mbr_lanczos_coeffs(mbr_lanczos *, double *, double *, void *) { MBR_FAIL(MBR_EUNSUPPORTED, "not built"); }
mbr_status mbr_lanczos_destroy(mbr_lanczos *) { return MBR_OK; }
mbr_status mbr_tridiag_lowest(const double *, const double *, const int32_t *, int32_t, int32_t, double *, void *) { MBR_FAIL(MBR_EUNSUPPORTED, "not built"); }
}
