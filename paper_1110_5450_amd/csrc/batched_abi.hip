// batched_abi.hip -- batched evaluation and the adjoint (C ABI).
#include <hip/hip_runtime.h>

#include "abi_internal.hpp"

using namespace sweep;

extern "C" {

size_t sweep_batched_workspace_size(const sweep_batch* batch, const sweep_options* opt) { (void)batch; (void)opt; return 0; }

sweep_status sweep_eval_batched(const sweep_batch* batch, const sweep_options* opt, void* pos, void* nrm,
                                void* workspace, size_t ws_bytes, void* stream)
{
    (void)batch; (void)opt; (void)pos; (void)nrm; (void)workspace; (void)ws_bytes; (void)stream;
    return fail(SWEEP_ERR_UNSUPPORTED, "not built yet");
}

size_t sweep_backward_workspace_size(const sweep_batch* batch, const sweep_options* opt) { (void)batch; (void)opt; return 0; }

sweep_status sweep_backward(const sweep_batch* batch, const sweep_options* opt, const void* grad_pos,
                            double* grad_path_ctrl, double* grad_prof_ctrl, void* workspace, size_t ws_bytes,
                            void* stream)
{
    (void)batch; (void)opt; (void)grad_pos; (void)grad_path_ctrl; (void)grad_prof_ctrl; (void)workspace; (void)ws_bytes; (void)stream;
    return fail(SWEEP_ERR_UNSUPPORTED, "not built yet");
}

void sweep_release_caches(void) {}

}
