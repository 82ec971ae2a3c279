// pending.hip -- entry points whose implementation lands in later files.
#include "../../include/mlspgemm.h"

extern "C" {

spgemm_status spgemm_batch_plan_create(int32_t, const spgemm_csr *, const spgemm_csr *, spgemm_csr *, int32_t, int32_t,
                                       void *, size_t, hipStream_t, spgemm_batch_plan **) { return SPGEMM_ERR_UNSUPPORTED; }
spgemm_status spgemm_batch_plan_run(spgemm_batch_plan *, hipStream_t) { return SPGEMM_ERR_UNSUPPORTED; }
void spgemm_batch_plan_destroy(spgemm_batch_plan *) {}

}
