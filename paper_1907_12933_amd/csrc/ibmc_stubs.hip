// Entry points whose kernels are not built yet report IBMC_E_UNIMPL.
#include "ibmc_host.h"

using namespace ibmc;

#define IBMC_STUB(name)                                                                           \
    return fail(IBMC_E_UNIMPL, #name " is not available in this build")

extern "C" ibmc_status ibmc_coverage(ibmc_ctx *, const ibmc_mlp *, const uint8_t *, const uint8_t *, int64_t, int32_t,
                                     const ibmc_cov_params *, ibmc_cov_summary *, uint64_t *) { IBMC_STUB(ibmc_coverage); }
extern "C" ibmc_status ibmc_coverage_dev(ibmc_ctx *, const ibmc_mlp *, const uint8_t *, const uint8_t *, int64_t,
                                         int32_t, const ibmc_cov_params *, ibmc_cov_summary *, uint64_t *) {
    IBMC_STUB(ibmc_coverage_dev);
}
extern "C" ibmc_status ibmc_coverage_all_dev(ibmc_ctx *, const ibmc_mlp *, const uint8_t *, const uint8_t *, int64_t,
                                             const ibmc_cov_params *, ibmc_cov_summary *, uint64_t *) {
    IBMC_STUB(ibmc_coverage_all_dev);
}
extern "C" ibmc_status ibmc_coverage_from_potentials(ibmc_ctx *, int32_t, const int32_t *, const int64_t *,
                                                     const int64_t *, int64_t, int32_t, const ibmc_cov_params *,
                                                     ibmc_cov_summary *, uint64_t *) {
    IBMC_STUB(ibmc_coverage_from_potentials);
}
extern "C" ibmc_status ibmc_proposer_create(ibmc_ctx *, uint64_t, ibmc_proposer **) { IBMC_STUB(ibmc_proposer_create); }
extern "C" void ibmc_proposer_free(ibmc_proposer *) {}
extern "C" ibmc_status ibmc_proposer_get(ibmc_proposer *, float *, float *, float *, float *) { IBMC_STUB(ibmc_proposer_get); }
extern "C" ibmc_status ibmc_proposer_set(ibmc_proposer *, const float *, const float *, const float *, const float *) {
    IBMC_STUB(ibmc_proposer_set);
}
extern "C" ibmc_status ibmc_proposer_features(ibmc_ctx *, const ibmc_mlp *, const uint8_t *, int32_t, int32_t,
                                              const int16_t *, int32_t, float *) { IBMC_STUB(ibmc_proposer_features); }
extern "C" ibmc_status ibmc_proposer_grad(ibmc_ctx *, ibmc_proposer *, const float *, const float *, int32_t, float,
                                          float *, float *, float *, float *, float *) { IBMC_STUB(ibmc_proposer_grad); }
extern "C" ibmc_status ibmc_proposer_train(ibmc_ctx *, ibmc_proposer *, const float *, const float *, int64_t,
                                           const ibmc_train_opts *, float *) { IBMC_STUB(ibmc_proposer_train); }
extern "C" ibmc_status ibmc_proposer_score(ibmc_ctx *, const ibmc_proposer *, const ibmc_mlp *, const uint8_t *,
                                           int32_t, int32_t, const int16_t *, int32_t, float *) {
    IBMC_STUB(ibmc_proposer_score);
}
extern "C" ibmc_status ibmc_check_property_ranked(ibmc_ctx *, const ibmc_mlp *, const ibmc_proposer *,
                                                  const uint8_t *, int32_t, int32_t, int32_t, const int16_t *, int32_t,
                                                  const ibmc_check_opts *, ibmc_check_summary *, ibmc_cex *) {
    IBMC_STUB(ibmc_check_property_ranked);
}
extern "C" ibmc_status ibmc_autotune(ibmc_ctx *, const ibmc_mlp *, int32_t, int32_t, char *, int64_t) {
    IBMC_STUB(ibmc_autotune);
}
