// Entry points that are not part of the plain forward path yet.
#include <hip/hip_runtime.h>

#include "dis.h"
#include "dis_host.h"

struct BatchPlan {
    int dummy;
};

void dis_batch_plan_free(BatchPlan* bp) { delete bp; }

extern "C" int dis_compute_flow_batched(dis_handle* h, int, const void* const*, const void* const*, const int*,
                                        const int*, const int*, void* const*) {
    if (!h) return DIS_EINVAL;
    h->err = "batched flow not built yet";
    return DIS_ESTATE;
}

extern "C" int dis_flow_backward(dis_handle* h, const void*, void*, void*) {
    if (!h) return DIS_EINVAL;
    h->err = "backward not built yet";
    return DIS_ESTATE;
}

extern "C" int dis_autotune(dis_handle* h, const char*) {
    if (!h) return DIS_EINVAL;
    return DIS_OK;
}
