// a5: batched form (placeholder until the persistent batched scheduler lands).
#include "common.h"

struct pardtw_plan {
    int32_t batch;
};

extern "C" pardtw_status pardtw_plan_create(int32_t batch, const int64_t* n_host, const int64_t* m_host, int64_t d,
                                            pardtw_prec prec, pardtw_plan** plan) {
    (void)batch; (void)n_host; (void)m_host; (void)d; (void)prec;
    if (plan) *plan = nullptr;
    return PARDTW_ERR_UNSUPPORTED;
}
extern "C" size_t pardtw_plan_workspace_bytes(const pardtw_plan* plan) { (void)plan; return 0; }
extern "C" int64_t pardtw_plan_path_capacity(const pardtw_plan* plan) { (void)plan; return 0; }
extern "C" void pardtw_plan_destroy(pardtw_plan* plan) { delete plan; }
extern "C" pardtw_status pardtw_align_batch(const pardtw_plan*, const float*, const float*, void*, size_t, float*,
                                            int32_t*, int32_t*, int32_t*, hipStream_t) {
    return PARDTW_ERR_UNSUPPORTED;
}
extern "C" pardtw_status pardtw_path_grad_batch(const pardtw_plan*, const float*, const float*, const int32_t*,
                                                const int32_t*, const float*, float*, float*, hipStream_t) {
    return PARDTW_ERR_UNSUPPORTED;
}
