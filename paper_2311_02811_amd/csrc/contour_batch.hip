// contour_batch.hip -- batched solve of many independent graphs.
#include <hip/hip_runtime.h>

#include "contour.h"
#include "contour_runtime.hpp"

extern "C" {

int contour_batch_plan_create(const contour_batch_t* batch, const contour_opts_t* opts,
                              contour_plan_t* plan_out)
{
    (void)batch;
    (void)opts;
    if (plan_out) *plan_out = nullptr;
    return CONTOUR_ENOTSUP;
}

int contour_batch_plan_launch(contour_plan_t plan, contour_stream_t stream)
{
    (void)plan;
    (void)stream;
    return CONTOUR_ENOTSUP;
}

int contour_batch_plan_destroy(contour_plan_t plan)
{
    (void)plan;
    return CONTOUR_OK;
}

int contour_cc_batched(const contour_batch_t* batch, const contour_opts_t* opts, contour_stream_t stream)
{
    (void)batch;
    (void)opts;
    (void)stream;
    return CONTOUR_ENOTSUP;
}

}  // extern "C"
