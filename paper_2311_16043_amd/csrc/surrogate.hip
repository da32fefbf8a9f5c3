// surrogate.hip -- MLP visibility surrogate (placeholder entry points).
#include "rv_internal.h"

using namespace rv;

extern "C" size_t rv_surrogate_bytes(void) { return 0; }
extern "C" size_t rv_surrogate_train_workspace_bytes(int32_t) { return 0; }
extern "C" size_t rv_surrogate_infer_workspace_bytes(int64_t) { return 0; }
extern "C" rv_status rv_surrogate_init(void *, uint64_t, const float *, const float *, void *) {
    set_error("rv_surrogate_init: not implemented");
    return RV_ERR_UNSUPPORTED;
}
extern "C" rv_status rv_surrogate_train(void *, const float *, const float *, const float *, int64_t,
                                        const rv_train_opts *, float *, void *, size_t, void *) {
    set_error("rv_surrogate_train: not implemented");
    return RV_ERR_UNSUPPORTED;
}
extern "C" rv_status rv_surrogate_infer_xd(const void *, const float *, const float *, int64_t, float *, float *,
                                           void *) {
    set_error("rv_surrogate_infer_xd: not implemented");
    return RV_ERR_UNSUPPORTED;
}
extern "C" rv_status rv_surrogate_infer(const void *, const void *, const rv_gaussians *, const float *, int32_t,
                                        const rv_trace_params *, int64_t, int64_t, float, float *, float *,
                                        int64_t *, void *, size_t, void *) {
    set_error("rv_surrogate_infer: not implemented");
    return RV_ERR_UNSUPPORTED;
}
