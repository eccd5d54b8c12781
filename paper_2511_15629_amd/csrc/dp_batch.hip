// Batched solves (placeholder until the persistent batched kernel lands).
#include "dpgpu.h"

struct dp_batch_plan {
    int n;
};

extern "C" {

int dp_batch_plan_create(dp_batch_plan **out, int n, const dp_problem *probs,
                         const char *tune_cache, void *stream)
{
    (void)out; (void)n; (void)probs; (void)tune_cache; (void)stream;
    return DP_ENOTSUP;
}

int dp_batch_solve(dp_batch_plan *plan, const float *const *lam, const float *const *P,
                   float *const *V1, int16_t *const *policy, void *stream)
{
    (void)plan; (void)lam; (void)P; (void)V1; (void)policy; (void)stream;
    return DP_ENOTSUP;
}

int dp_batch_solve_looped(dp_batch_plan *plan, const float *const *lam, const float *const *P,
                          float *const *V1, int16_t *const *policy, void *stream)
{
    (void)plan; (void)lam; (void)P; (void)V1; (void)policy; (void)stream;
    return DP_ENOTSUP;
}

int dp_batch_plan_describe(const dp_batch_plan *plan, char *buf, size_t len)
{
    (void)plan; (void)buf; (void)len;
    return DP_ENOTSUP;
}

void dp_batch_plan_destroy(dp_batch_plan *plan) { (void)plan; }

}
