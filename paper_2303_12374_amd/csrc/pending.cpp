// Batched and served forms: entry points present, implementation pending.
#include "kl_internal.hpp"

using namespace kl;

extern "C" {
int kl_batch_create(const kl_grid_t *, void *const *, int32_t, double, int32_t, void *, void **)
{
    return fail(KL_ERR_INVALID, "batched form not available in this build");
}
int kl_batch_run(void *, void *) { return fail(KL_ERR_INVALID, "batched form not available"); }
int kl_batch_info(void *, int32_t *, int64_t *) { return fail(KL_ERR_INVALID, "batched form not available"); }
int kl_batch_destroy(void *) { return fail(KL_ERR_INVALID, "batched form not available"); }
int kl_server_create(void *, size_t, size_t, void **) { return fail(KL_ERR_INVALID, "server not available"); }
int kl_submit(void *, const kl_request_t *, uint64_t *) { return fail(KL_ERR_INVALID, "server not available"); }
int kl_poll(void *, uint64_t, kl_result_t *) { return fail(KL_ERR_INVALID, "server not available"); }
int kl_release(void *, uint64_t) { return fail(KL_ERR_INVALID, "server not available"); }
int kl_server_stats(void *, int64_t *) { return fail(KL_ERR_INVALID, "server not available"); }
int kl_server_destroy(void *) { return fail(KL_ERR_INVALID, "server not available"); }
}
