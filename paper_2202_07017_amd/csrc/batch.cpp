// Batched evaluation of many small rotation circuits (energies and adjoint
// gradients) -- placeholder entry points until the persistent kernel lands.
#include "qsv.h"
#include "qsv_host.h"

using namespace qsv;

struct qsv_batch_plan {
    int ninst = 0;
};

extern "C" {

qsv_status qsv_batch_plan_create(const qsv_circuit*, const qsv_pauli_sum*, int, qsv_dtype,
                                 qsv_batch_plan**, size_t*)
{
    return fail(QSV_ERR_UNSUPPORTED, "batched evaluation is not available in this build");
}

qsv_status qsv_batch_offsets(const qsv_batch_plan*, int64_t*)
{
    return fail(QSV_ERR_UNSUPPORTED, "batched evaluation is not available in this build");
}

qsv_status qsv_batch_run(qsv_batch_plan*, const double*, void*, double*, double*, void*)
{
    return fail(QSV_ERR_UNSUPPORTED, "batched evaluation is not available in this build");
}

qsv_status qsv_batch_tune(qsv_batch_plan*, const double*, void*, double*, double*, void*, int*)
{
    return fail(QSV_ERR_UNSUPPORTED, "batched evaluation is not available in this build");
}

qsv_status qsv_batch_plan_destroy(qsv_batch_plan* plan)
{
    delete plan;
    return ok();
}

}  // extern "C"
