// grad.hip -- reverse mode of the deterministic stream (see psvd.h).
#include <hip/hip_runtime.h>

#include "kernels.h"

extern "C" int psvd_stream_backward(const void*, int64_t, int64_t, int32_t, int32_t, int64_t, int32_t, double,
                                    const void*, const double*, void*, void*) {
    return PSVD_E_STATE;
}

extern "C" int psvd_loss_grad(const void*, int64_t, int64_t, int32_t, int32_t, int64_t, int32_t, double,
                              const double*, double*, void*, void*) {
    return PSVD_E_STATE;
}
